"""CPU FP64 oracle for non-zero noise extrapolation (arxiv 2501.13237).

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
executes anything in this directory; only ``tests/``, the smoke check in
``__graft_entry__.py`` and the ``cpu_baseline`` leg of ``bench.py`` use it.

The oracle is a plain, slow, obviously correct restatement of what the paper's
method computes, written in NumPy float64 / complex128:

* ``ptm``       -- Pauli-transfer matrices of gates and noise channels
                   (Sec. 2.2.1 "Parametrised noise models", App. C.2).
* ``dense``     -- brute-force 2^n x 2^n density-matrix simulation with Kraus
                   operators in the computational basis (independent check).
* ``pauliprop`` -- exact Heisenberg-picture Pauli propagation for Clifford
                   gates under Pauli noise (independent check).
* ``mpo``       -- the vectorised-MPO emulation of Sec. 2.1 in the real Pauli
                   basis: zig-zag two-site updates, truncated SVD to a fixed
                   bond dimension, partial/emulation fidelity, readout.
* ``mpo_ketbra``-- the same emulation in the paper's complex ket-bra superket
                   basis (eq. ``vectorized_dm``), used to pin the Pauli-basis
                   oracle by basis invariance.
* ``fits``      -- the noise-strength extrapolations of Sec. 2.2.2 (B) and
                   App. B.2, the polynomial fit, and the fidelity
                   extrapolation of Sec. 2.2.2 (A) with App. B.1's criterion.

It shares no code with the HIP/C++ path.
"""
