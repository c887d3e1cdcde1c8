"""The tuner: it measures launch parameters on the device and MPOs created
with block = 0 follow its record.  Group size and kernel build never change a
result (bitwise); the cross-block-only schedule changes the rotation order,
so those results agree with the defaults within the path's tolerance."""
import sys

import numpy as np
import pytest

from oracle import mpo as ompo
from oracle import ptm
from paper_2501_13237_amd import nze, workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(n, chi, layers, noise, factors, precision, block):
    m = nze.MPO(n, chi, len(factors), precision, block=block)
    nze.run_circuit(m, layers, noise, factors)
    out = m.expect(workloads.z_singles(n) + workloads.zz_neighbours(n))
    m.close()
    return out


@pytest.mark.parametrize("precision,tol", [(nze.NZE_FP64, 1e-10), (nze.NZE_MIXED, 1e-5)])
def test_tuned_launches_match_defaults(precision, tol):
    n, chi = 14, 64
    factors = [1.0, 2.0, 4.0, 8.0]
    noise = {"dep": 2e-3}
    layers = workloads.brickwork(n, 10, seed=71)
    rec = nze.tune(chi, precision, len(factors))
    _say(f"tuned prec={precision}: {rec}")
    assert rec["block"] == 16 and rec["group_scale"] in (1, 2) and rec["kernel"] in (1, 2)
    assert rec["ms_per_svd"] > 0 and nze.tuning_get(chi, precision, len(factors)) == rec
    ref = _run(n, chi, layers, noise, factors, precision, 16)
    got = _run(n, chi, layers, noise, factors, precision, 0)
    if (rec["cross_sweeps"], rec["cross_min_blocks"]) == (8, 64):
        assert all(np.array_equal(a, b) for a, b in zip(ref, got))
    # every launch choice with the default schedule is bitwise the default
    for scale in (1, 2):
        for kernel in ((1, 2) if precision == nze.NZE_MIXED else (1,)):
            nze.tuning_set(chi, precision, len(factors),
                           dict(block=16, group_scale=scale, kernel=kernel, cross_sweeps=8,
                                cross_min_blocks=64, ms_per_svd=1.0))
            got = _run(n, chi, layers, noise, factors, precision, 0)
            assert all(np.array_equal(a, b) for a, b in zip(ref, got)), (scale, kernel)
    # another schedule: within tolerance of the defaults and of the oracle
    nze.tuning_set(chi, precision, len(factors),
                   dict(block=16, group_scale=1, kernel=1, cross_sweeps=4,
                        cross_min_blocks=16, ms_per_svd=1.0))
    got = _run(n, chi, layers, noise, factors, precision, 0)
    assert np.max(np.abs(got[0] - ref[0])) < tol
    obs = workloads.z_singles(n) + workloads.zz_neighbours(n)
    for j, c in enumerate(factors):
        m = ompo.PauliMPO(n, chi, tie_tol=1e-10 if precision == nze.NZE_FP64 else 1e-5)
        nz = ptm.Noise(**noise).scaled(c)
        for ls, us in layers:
            m.apply_layer(ls, [ptm.ptm_noisy_gate(U, nz) for U in us])
        assert np.max(np.abs(got[0][j] - m.expectations(obs))) < tol
    nze.tuning_set(chi, precision, len(factors), rec)
