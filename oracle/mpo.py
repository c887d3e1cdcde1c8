"""Vectorised-MPO emulation of a noisy circuit in the real Pauli basis.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

What is computed (paper Sec. 2.1):

* State representation (Sec. 2.1.1): the vectorised density operator is an MPS
  of local dimension 4 and bond dimension at most D (here ``chi_max``).  Site k
  holds M[k] of shape (chi_left, 4, chi_right).  The local index is the Pauli
  coordinate v_P = Tr(P rho) (P in I, X, Y, Z), a fixed orthogonal change of
  basis (up to a factor sqrt(2) per site) of the paper's ket-bra superket index
  (i_k, j_k), so singular values, truncations, fidelities and expectation
  values are the same in both bases (pinned by ``oracle.mpo_ketbra``).
* Approximate emulation (Sec. 2.1.2): one subcircuit C_l is one noisy
  two-qubit gate.  C_l is applied to the current approximate state and the
  result is replaced by the closest (Frobenius) state of bond dimension at most
  D, renormalised to Frobenius norm 1; the initial state is a product state.
  The closest state is obtained, as usual, by bringing the MPO into mixed
  canonical form around the two sites of the gate (App. A.1's footnote on
  canonical form), contracting the two sites, applying the gate's 16x16
  superoperator and truncating the SVD of the two-site block.
* Partial fidelity (Sec. 2.1.2, eq. for f_l): with orthonormal environments the
  two-site block carries the whole state, the truncation is the orthogonal
  projection onto the leading singular vectors, and f_l reduces to
  (sum of kept s_i^2) / (sum of all s_i^2).  The emulation fidelity is the
  product of the f_l (eq. ``emulation_fidelity``).
* Readout: <P> = Tr(P rho) / Tr(rho) = c_P / c_I, where c_X is the contraction
  of the Pauli-X_k slices of every site ("up to normalization", Sec. 2.1.2).

Readings where the paper is silent (recorded in the design notes):

* Schedule: the gates of one layer are applied one at a time in zig-zag
  order -- increasing left site when the layer's left sites are even (left to
  right), decreasing when they are odd (right to left).  Before a gate on
  (k, k+1) the orthogonality centre is moved to k (left to right) or k+1
  (right to left) by QR / LQ steps.  After a left-to-right gate the new M[k] is
  U_r (left-orthonormal) and M[k+1] = S_r V_r^T; right to left, M[k] = U_r S_r
  and M[k+1] = V_r^T.
* Truncation rule: r = min(chi_max, #{s_i > tau * s_1}), r >= 1.  If the cut is
  set by chi_max and the last kept and first dropped values agree within
  relative ``tie_tol``, the whole (chained) cluster of tied values is dropped;
  if that would drop everything, r = chi_max.
* Normalisation: the centre is renormalised to Frobenius norm 1 after every
  gate and the logarithm of the removed factor is accumulated in
  ``log_scale``, so exp(log_scale) * c_I is the trace of the (truncated) state.
"""
import numpy as np


def truncation_rank(s, chi_max, tau, tie_tol):
    """Number of singular values kept (``s`` sorted in decreasing order)."""
    s = np.asarray(s, dtype=np.float64)
    if s.size == 0 or s[0] <= 0.0:
        return 1
    above = int(np.count_nonzero(s > tau * s[0]))
    r = max(1, min(chi_max, above))
    if r == chi_max and r < above:
        r0 = r
        while r > 0 and (s[r - 1] - s[r]) <= tie_tol * s[r - 1]:
            r -= 1
        if r == 0:
            r = r0
    return r


def product_site(bit):
    """Pauli coordinates (Tr(I rho), Tr(X rho), Tr(Y rho), Tr(Z rho)) of
    |bit><bit|."""
    return np.array([1.0, 0.0, 0.0, -1.0 if bit else 1.0])


class PauliMPO:
    def __init__(self, n, chi_max, tau=1e-14, tie_tol=1e-10, init_bits=None,
                 init_sites=None):
        self.n = n
        self.chi_max = chi_max
        self.tau = tau
        self.tie_tol = tie_tol
        if init_sites is None:
            bits = init_bits if init_bits is not None else [0] * n
            init_sites = [product_site(b) for b in bits]
        self.sites = []
        self.log_scale = 0.0
        for v in init_sites:
            v = np.asarray(v, dtype=np.float64)
            nv = np.linalg.norm(v)
            self.sites.append((v / nv).reshape(1, 4, 1))
            self.log_scale += np.log(nv)
        self.centre = 0
        self.fidelity = 1.0
        self.partial_fidelities = []
        self.discarded = []          # discarded weight 1 - f per gate
        self.cut_gaps = []           # relative gap (s_r - s_{r+1}) / s_1 at cuts

    # ------------------------------------------------------------ canonical
    def move_centre(self, target):
        """QR (left to right) / LQ (right to left) steps, one site at a time."""
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
            Q, R = np.linalg.qr(M.reshape(cl, 4 * cr).T)   # M = R^T Q^T
            self.sites[c] = Q.T.reshape(Q.shape[1], 4, cr)
            self.sites[c - 1] = np.einsum('apj,jk->apk', self.sites[c - 1],
                                          R.T)
            self.centre -= 1

    # ------------------------------------------------------------- updates
    def two_site_block(self, k, R):
        """Theta' = (R x 1) Theta as a (4 chi_l) x (4 chi_r) matrix, rows
        (a, p'), columns (q', b)."""
        A, B = self.sites[k], self.sites[k + 1]
        cl, cr = A.shape[0], B.shape[2]
        theta = np.einsum('apc,cqb->apqb', A, B).reshape(cl, 16, cr)
        theta = np.einsum('PQ,aQb->aPb', R, theta)
        return theta.reshape(cl * 4, 4 * cr)

    def apply_gate(self, k, R, left_to_right):
        self.move_centre(k if left_to_right else k + 1)
        cl, cr = self.sites[k].shape[0], self.sites[k + 1].shape[2]
        Xm = self.two_site_block(k, np.asarray(R, dtype=np.float64))
        try:
            U, s, Vt = np.linalg.svd(Xm, full_matrices=False)
        except np.linalg.LinAlgError:
            import scipy.linalg
            U, s, Vt = scipy.linalg.svd(Xm, full_matrices=False,
                                        lapack_driver='gesvd')
        r = truncation_rank(s, self.chi_max, self.tau, self.tie_tol)
        s2 = s * s
        kept, total = s2[:r].sum(), s2.sum()
        f = kept / total
        if r < s.size:
            self.cut_gaps.append((s[r - 1] - s[r]) / s[0])
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
        self.discarded.append(1.0 - f)
        return f

    def apply_layer(self, left_sites, ptms):
        """Apply one layer of gates on pairs (k, k+1), k in ``left_sites``
        (strictly increasing, pairs disjoint), ``ptms[i]`` being the 16x16
        superoperator of the gate on ``left_sites[i]``."""
        ls = list(left_sites)
        if any(b - a < 2 for a, b in zip(ls, ls[1:])):
            raise ValueError("left sites must be increasing and disjoint")
        if ls and (ls[0] < 0 or ls[-1] + 1 >= self.n):
            raise ValueError("gate outside the chain")
        if not ls:
            return
        ltr = (ls[0] % 2 == 0)
        order = range(len(ls)) if ltr else range(len(ls) - 1, -1, -1)
        for i in order:
            self.apply_gate(ls[i], ptms[i], ltr)

    # ------------------------------------------------------------- readout
    def contract(self, paulis):
        v = np.ones(1)
        for k, p in enumerate(paulis):
            v = v @ self.sites[k][:, int(p), :]
        return v[0]

    def expectations(self, observables):
        cI = self.contract([0] * self.n)
        return np.array([self.contract(o) / cI for o in observables])

    def trace(self):
        return np.exp(self.log_scale) * self.contract([0] * self.n)

    def bond_dims(self):
        return [self.sites[k].shape[2] for k in range(self.n - 1)]

    def bond_spectrum(self, l):
        """Schmidt values across bond (l, l+1) of the normalised state."""
        saved = ([s.copy() for s in self.sites], self.centre)
        self.move_centre(l)
        M = self.sites[l]
        s = np.linalg.svd(M.reshape(M.shape[0] * 4, M.shape[2]),
                          compute_uv=False)
        self.sites, self.centre = saved
        return s

    def entanglement_entropy(self, l):
        """MPO entanglement entropy at bond l (App. A.1)."""
        s = self.bond_spectrum(l)
        p = s * s / np.sum(s * s)
        p = p[p > 0]
        return float(-np.sum(p * np.log(p)))

    def pauli_vector(self):
        """Full 4^n Pauli-coordinate vector v_P = Tr(P rho) (small n only)."""
        v = np.ones((1, 1))
        for M in self.sites:
            v = np.einsum('xa,apb->xpb', v, M).reshape(-1, M.shape[2])
        return np.exp(self.log_scale) * v[:, 0]


def run(n, layers, chi_max, tau=1e-14, tie_tol=1e-10, init_bits=None):
    """Evolve the product state through ``layers``, a list of
    (left_sites, ptms) pairs."""
    m = PauliMPO(n, chi_max, tau, tie_tol, init_bits=init_bits)
    for left_sites, ptms in layers:
        m.apply_layer(left_sites, ptms)
    return m
