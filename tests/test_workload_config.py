"""The committed workload configuration (synth/workloads.json) is the
module's, and its method constants are the ones the code uses."""
import inspect
import json
import math
import os

from synth import cluster as SC
from synth import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_json_matches_module():
    with open(os.path.join(ROOT, "synth", "workloads.json")) as f:
        assert json.load(f) == json.loads(json.dumps(W.as_config()))


def test_method_constants_match_the_code():
    m = W.METHOD
    from paper_2303_00790_amd import scf
    d = {k: v.default for k, v in inspect.signature(scf.setup).parameters.items()}
    assert d["margin"] == m["domain_margin_bohr"]
    assert d["mix_beta"] == m["anderson_beta"] and d["mix_history"] == m["anderson_history"]
    assert d["first_iters"] == m["chfsi_iters_first_scf_step"]
    assert SC.D_SIH == m["bond_si_h_angstrom"]
    assert SC.A_SI_OBSERVED == m["lattice_angstrom"] and SC.A_SI_OPTIMISED == m["lattice_table_i_angstrom"]
    for ne in (8, 142, 4121 * 2, 7000):
        assert SC.n_states(ne) == 64 * math.ceil(math.ceil(1.1 * ne / 2) / 64)
