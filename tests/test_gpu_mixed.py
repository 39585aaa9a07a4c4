"""Mixed precision: the FP32 filter (H X recurrences) and FP32-input MFMA Gram
products with FP64 Cholesky, eigensolve and mixing, run to self-consistency
and compared with the FP64 path (itself parity-tested against the oracle to
1e-8 Ha) from the same seed.  Bounds: 1e-5 Ha on the occupied eigenvalues and
1e-5 Ha per atom on the total energy."""
import numpy as np
import pytest

from synth.cluster import make_cluster
from synth.workloads import MODEL_PP

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _converge(dtype):
    from paper_2303_00790_amd import scf as S
    c = make_cluster(5.5, 1001)
    st = S.setup(c, MODEL_PP, dtype=dtype)
    rho0 = st["H"].sad_density(c.pos, c.species, c.n_electrons)
    res = S.run(st, rho0, max_steps=40, sre_tol_ry=1e-5)
    return c, res


def test_mixed_precision_matches_fp64():
    c, r64 = _converge("f64")
    _, r32 = _converge("f32")
    assert r64.converged and r32.converged, (r64.steps, r32.steps)
    occ = c.n_electrons // 2
    d_eig = np.abs(r32.eig[:occ] - r64.eig[:occ]).max()
    d_e = abs(r32.energy - r64.energy) / c.n_atoms
    print(f"mixed vs FP64: max |d eig| = {d_eig:.2e} Ha, |dE|/atom = {d_e:.2e} Ha, steps {r32.steps} vs {r64.steps}")
    assert d_eig < 1e-5
    assert d_e < 1e-5
    assert r64.reports[-1]["lumo"] - r64.reports[-1]["homo"] > 0.05
