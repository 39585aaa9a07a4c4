"""The trained initial-density network against the plain superposition start,
through the C ABI: both FP64 SCFs (same start vectors, the paper's schedule
of four ChFSI iterations then one, SRE < 1e-4 Ry) on one cluster the network
never saw (the record's test cluster: 2.5 nm, a geometry seed outside the
training seeds), the learned start from the committed weights (32-channel
network, its correction high-passed at 8 cells).

The learned start must take fewer SCF steps and reach the same energy within
1e-5 Ha per atom (the mixed-precision energy bound; both runs here are FP64,
so their converged energies differ only by where each stops).
"""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "results", "dnet_c32.npy")
RECORD = os.path.join(ROOT, "results", "learned_density_4nm.json")


def test_learned_start_saves_scf_steps():
    from paper_2303_00790_amd import binding as B
    from paper_2303_00790_amd import density_model as DM
    from synth.cluster import make_cluster
    from synth.workloads import MODEL_PP
    rec = json.load(open(RECORD))
    case = rec["test_cluster"]
    net = B.DensityNet(rec["channels"], seed=1)
    net.set_params(np.load(WEIGHTS).astype(np.float32))
    c = make_cluster(5.0 * case["diam_nm"], case["seed"], sigma_angstrom=0.02)
    row = DM.evaluate(net, [c], MODEL_PP, dtype="f64", highpass_sigma=rec["highpass_sigma"],
                      log=lambda m: print(m, flush=True))[0]
    print(row)
    assert row["conv_sad"] and row["conv_net"]
    assert row["steps_net"] < row["steps_sad"], row
    assert row["de_per_atom"] <= 1e-5, row
