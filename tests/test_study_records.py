"""Host logic of the study drivers (CPU): the mixed-vs-FP64 comparison
record, the merge of density-network training and evaluation records, and
the merge and refit of gap-study runs, on hand-made records whose results
are known."""
import json

import numpy as np
import pytest

from paper_2303_00790_amd import gap_study, precision_study, train_density


def test_precision_compare_reports_differences_of_the_two_runs():
    info = dict(workload="w", n_si=3, n_h=1, n_atoms=4, degree=12)
    r64 = dict(eig_occ=[-1.0, -0.5, -0.25], energy=-10.0, steps=10, seconds=20.0, n_points=100, M=64,
               sre_tol=1e-5, sre_last=5e-6, converged=True, start_density="rho.npy")
    r32 = dict(eig_occ=[-1.0 + 2e-6, -0.5 - 4e-6, -0.25], energy=-10.0 + 8e-6, steps=8, seconds=8.0,
               n_points=100, M=64, sre_tol=1e-5, sre_last=7e-6, converged=True, start_density="rho.npy")
    c = precision_study.compare(info, r64, r32)
    assert c["max_occ_eig_diff_ha"] == pytest.approx(4e-6)
    assert c["mean_occ_eig_diff_ha"] == pytest.approx(2e-6)
    assert c["de_per_atom_ha"] == pytest.approx(2e-6)
    assert c["s_per_step_f64"] == 2.0 and c["s_per_step_mixed"] == 1.0
    assert c["start_density_f64"] == c["start_density_mixed"] == "rho.npy"
    assert c["converged"]
    r32["converged"] = False
    assert not precision_study.compare(info, r64, r32)["converged"]


def _eval(seeds, steps, diam=4.0):
    rows = [dict(n_atoms=100, steps_sad=a, steps_net=b, conv_sad=True, conv_net=True, e_sad=-1.0, e_net=-1.0,
                 de_per_atom=1e-9 * (i + 1), sre0_sad=10.0, sre0_net=5.0) for i, (a, b) in enumerate(steps)]
    return dict(channels=32, dtype="f64", eval_diam_nm=diam, eval_seeds=seeds, first_iters=4, highpass_sigma=8.0,
                eval=rows)


def test_density_records_merge(tmp_path):
    train = dict(channels=32, dtype="f64", train_clusters=120, steps=2000, patch=64, loss_first=0.3, loss_last=0.01)
    paths = []
    for name, rec in (("t", train), ("a", _eval([1, 2], [(40, 30), (38, 34)])), ("b", _eval([3], [(42, 32)]))):
        p = tmp_path / f"{name}.json"
        p.write_text(json.dumps(rec))
        paths.append(str(p))
    tp = tmp_path / "test.json"
    tp.write_text(json.dumps(_eval([9], [(25, 21)], diam=2.5)))
    res = train_density.merge_records(paths, str(tp))
    assert res["eval_seeds"] == [1, 2, 3]
    assert res["mean_steps_sad"] == pytest.approx(40.0)
    assert res["mean_steps_net"] == pytest.approx(32.0)
    assert res["max_de_per_atom"] == pytest.approx(2e-9)
    assert res["train"]["train_clusters"] == 120
    assert res["test_cluster"] == dict(diam_nm=2.5, seed=9, highpass_sigma=8.0, dtype="f64", steps_sad=25,
                                       steps_net=21, de_per_atom=1e-9)
    assert res["small_clusters"]["seeds"] == [9] and len(res["small_clusters"]["eval"]) == 1
    other = tmp_path / "c.json"
    other.write_text(json.dumps(_eval([4], [(40, 30)], diam=3.0)))
    with pytest.raises(SystemExit):
        train_density.merge_records(paths + [str(other)])


def test_gap_study_merge_refits_the_joined_clusters(tmp_path):
    # gaps on the curve E0 + A / d^k exactly: the free fit returns it
    e0, a, k = 1.1, 2.3, 1.4
    pp = dict(r_loc=0.7)
    runs = []
    for ds in ((1.0, 2.0, 3.0), (4.0, 5.0)):
        rows = [dict(diam_nm=d, gap_ev=e0 + a / d ** k) for d in ds]
        p = tmp_path / f"g{len(runs)}.json"
        p.write_text(json.dumps(dict(h=0.7, dtype="f32", pp=pp, clusters=rows)))
        runs.append(str(p))
    out = tmp_path / "all.json"
    res = gap_study.main(["--merge", runs[1], runs[0], "--out", str(out)])
    assert [c["diam_nm"] for c in res["clusters"]] == [1.0, 2.0, 3.0, 4.0, 5.0]
    saved = json.loads(out.read_text())
    assert saved["fit"]["e0_ev"] == pytest.approx(e0, rel=1e-4)
    assert saved["fit"]["a_ev"] == pytest.approx(a, rel=1e-4)
    assert saved["fit"]["k"] == pytest.approx(k, rel=1e-4)
    bad = tmp_path / "bad.json"
    bad.write_text(json.dumps(dict(h=0.9, dtype="f32", pp=pp, clusters=[])))
    with pytest.raises(SystemExit):
        gap_study.main(["--merge", runs[0], str(bad)])
