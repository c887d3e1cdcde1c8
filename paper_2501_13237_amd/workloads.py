"""Seeded synthetic inputs: brickwork circuits, noise levels, observables.

This module generates inputs only and holds none of the method's arithmetic:
it produces 4x4 gate unitaries, noise parameters, amplification factors and
Pauli strings.  Both the library (through its C-ABI) and the test oracle take
these as inputs; neither builds them itself.

* Haar-random SU(4): QR of a complex Ginibre matrix with the phases of R's
  diagonal moved into Q (Mezzadri, "How to generate random matrices from the
  classical compact groups", 2007), then the determinant phase removed.
* Random two-qubit Clifford: uniform over the 11520 elements of the two-qubit
  Clifford group modulo global phase, enumerated once by breadth-first search
  from {H x I, I x H, S x I, I x S, CNOT}.
* Brickwork on a 1D open chain: layer t acts on pairs (k, k+1) with
  k = t (mod 2).
"""
from dataclasses import dataclass, field

import numpy as np

# ------------------------------------------------------------------ gates


def haar_su4(rng):
    z = (rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))
    z /= np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    q = q * (d / np.abs(d))[None, :]
    q /= np.linalg.det(q) ** 0.25
    return q


_CLIFFORDS = None


def _phase_key(U):
    flat = U.reshape(-1)
    i = int(np.argmax(np.abs(flat) > 1e-6))
    ph = flat[i] / abs(flat[i])
    V = U / ph
    key = np.rint(np.concatenate([V.real, V.imag]).reshape(-1) * 1e6)
    return key.astype(np.int64).tobytes(), V


def clifford_group2():
    """All 11520 two-qubit Cliffords modulo phase, as 4x4 unitaries, in a
    deterministic order."""
    global _CLIFFORDS
    if _CLIFFORDS is not None:
        return _CLIFFORDS
    H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
    S = np.array([[1, 0], [0, 1j]], dtype=np.complex128)
    I = np.eye(2, dtype=np.complex128)
    CX = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]],
                  dtype=np.complex128)
    gens = [np.kron(H, I), np.kron(I, H), np.kron(S, I), np.kron(I, S), CX]
    k0, e = _phase_key(np.eye(4, dtype=np.complex128))
    seen = {k0: e}
    order = [e]
    frontier = [e]
    while frontier:
        nxt = []
        for U in frontier:
            for g in gens:
                k, V = _phase_key(g @ U)
                if k not in seen:
                    seen[k] = V
                    order.append(V)
                    nxt.append(V)
        frontier = nxt
    _CLIFFORDS = order
    return order


def random_clifford2(rng):
    group = clifford_group2()
    return group[int(rng.integers(len(group)))]


# --------------------------------------------------------------- circuits


def brickwork_left_sites(n, t):
    return list(range(t % 2, n - 1, 2))


def brickwork(n, depth, seed, kind="haar"):
    """List of layers; each layer is (left_sites, [U per gate])."""
    rng = np.random.default_rng(seed)
    draw = haar_su4 if kind == "haar" else random_clifford2
    layers = []
    for t in range(depth):
        ls = brickwork_left_sites(n, t)
        layers.append((ls, [draw(rng) for _ in ls]))
    return layers


def n_gates(layers):
    return sum(len(ls) for ls, _ in layers)


# ------------------------------------------------------------ observables


def pauli_string(n, ops):
    """ops: dict site -> 'X'|'Y'|'Z' (or 1..3); returns uint8[n]."""
    code = {"I": 0, "X": 1, "Y": 2, "Z": 3}
    s = np.zeros(n, dtype=np.uint8)
    for k, p in ops.items():
        s[k] = code[p] if isinstance(p, str) else int(p)
    return s


def z_singles(n):
    return [pauli_string(n, {i: "Z"}) for i in range(n)]


def zz_neighbours(n):
    return [pauli_string(n, {i: "Z", i + 1: "Z"}) for i in range(n - 1)]


def weight1_all(n):
    return [pauli_string(n, {i: p}) for i in range(n) for p in "XYZ"]


def weight2_neighbours(n):
    return [pauli_string(n, {i: p, i + 1: q}) for i in range(n - 1)
            for p in "XYZ" for q in "XYZ"]


# -------------------------------------------------------------- workloads


@dataclass
class Workload:
    name: str
    n: int
    depth: int
    kind: str                      # "haar" | "clifford"
    noise: dict                    # base noise parameters (p0 etc.)
    factors: list                  # amplification factors c_j
    chi: int
    observables: list = field(default_factory=list)
    seed: int = 0

    def circuit(self):
        return brickwork(self.n, self.depth, self.seed, self.kind)


def plain_fp64_n8(seed=0):
    """n = 8 chain, depth-8 Haar SU(4) brickwork, two-qubit depolarizing
    p = 1e-3 amplified by {1, 2, 4, 8}, chi = 256 (exact at n = 8)."""
    n = 8
    return Workload("haar-n8-d8-dep1e-3-L4-chi256", n, 8, "haar",
                    {"dep": 1e-3}, [1.0, 2.0, 4.0, 8.0], 256,
                    z_singles(n) + zz_neighbours(n), seed)


def mixed_n32(chi=64, seed=0):
    """n = 32 chain, depth 20, depolarizing 1e-3 plus amplitude damping
    gamma = 5e-4 on each qubit, one noise level; all <Z_i>."""
    n = 32
    return Workload(f"haar-n32-d20-dep1e-3-ad5e-4-chi{chi}", n, 20, "haar",
                    {"dep": 1e-3, "ad": 5e-4}, [1.0], chi, z_singles(n), seed)


def noise_sweep_n50(seed=0, levels=8):
    """n = 50 chain, depth 24, 8 levels lambda_j = (1 + 15 j / 7) p0 with
    p0 = 1e-3, chi = 256; <Z_25> and <X_1 X_2>."""
    n = 50
    factors = [1.0 + 15.0 * j / (levels - 1) for j in range(levels)]
    obs = [pauli_string(n, {25: "Z"}), pauli_string(n, {1: "X", 2: "X"})]
    return Workload("haar-n50-d24-dep1e-3-L8-chi256", n, 24, "haar",
                    {"dep": 1e-3}, factors, 256, obs, seed)


def clifford_n64(seed=0):
    """n = 64 chain, depth 30 random two-qubit Cliffords, Pauli noise
    px = py = pz = 3e-4 on each qubit, factors {1, 4, 7, 10, 13, 16},
    chi = 512; all weight-1 and nearest-neighbour weight-2 Paulis."""
    n = 64
    return Workload("clifford-n64-d30-pauli3e-4-L6-chi512", n, 30, "clifford",
                    {"px": 3e-4, "py": 3e-4, "pz": 3e-4},
                    [1.0, 4.0, 7.0, 10.0, 13.0, 16.0], 512,
                    weight1_all(n) + weight2_neighbours(n), seed)
