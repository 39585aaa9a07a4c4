"""Cross-checks of the hand-transcribed fixtures in tests/golden against the
figures the paper derives from them in its text (Results section), so that a
slip in transcribing Table I fails here rather than inside another pin."""
from golden import table_i, text_figures

FIG = text_figures()
ROWS = table_i()


def test_six_rows_in_size_order():
    assert len(ROWS) == 6
    assert [r.diameter_nm for r in ROWS] == sorted(r.diameter_nm for r in ROWS)
    assert [r.n_si for r in ROWS] == sorted(r.n_si for r in ROWS)


def test_names_match_counts():
    for r in ROWS:
        assert r.name == f"Si{r.n_si}H{r.n_h}"


def test_largest_degrees_of_freedom():
    # grid points times states of the largest cluster, as the text states it (two digits)
    big = ROWS[-1]
    assert round(big.grid_points * big.states / 1e12, 1) == FIG["degrees_of_freedom_largest"] / 1e12


def test_largest_computed_fraction():
    big = ROWS[-1]
    assert round(100 * big.states / big.grid_points, 2) == FIG["computed_fraction_percent"]


def test_spacing_ratio_and_spacings():
    assert round((0.7 / 0.9) ** 3, 2) == FIG["spacing_size_ratio"]
    # the two largest clusters use h = 0.9 bohr, the rest h = 0.7 bohr
    assert [r.h_bohr for r in ROWS] == [0.7] * 4 + [0.9] * 2


def test_lattice_constants_within_one_percent():
    opt, obs = FIG["lattice_optimised_angstrom"], FIG["lattice_observed_angstrom"]
    assert abs(opt - obs) / obs < 0.01


def test_grid_points_fill_a_sphere_larger_than_the_cluster():
    # every domain holds the cluster: (4/3) pi (d/2)^3 / h^3 is below the printed count
    bohr_nm = 0.0529177
    for r in ROWS:
        cluster_points = 4.0 / 3.0 * 3.141592653589793 * (r.diameter_nm / 2 / bohr_nm) ** 3 / r.h_bohr ** 3
        assert cluster_points < r.grid_points < 3 * cluster_points


def test_gap_fit_constants_are_physical():
    # a positive offset below silicon's LDA-scale gap, and an exponent between the earlier
    # small-cluster fits (1.1 to 1.39) and the effective-mass limit of 2, as the text argues
    assert 0 < FIG["gap_offset_ev"] < 1.2 and 1.39 < FIG["gap_exponent"] < 2.0
    assert 0.99 < FIG["gap_fit_r2"] < 1.0


def test_oracle_scf_reference_is_consistent():
    # the computed fixture: occupied eigenvalues ascending, HOMO the last of
    # them, a gap to the LUMO, one state per electron pair, converged below
    # the threshold the generator uses
    import json
    from pathlib import Path
    ref = json.loads((Path(__file__).resolve().parent / "golden" / "scf_si35_oracle.json").read_text())
    e = ref["eig_occ_ha"]
    assert len(e) == ref["cluster"]["n_electrons"] // 2
    assert all(a <= b for a, b in zip(e, e[1:]))
    assert e[-1] == ref["homo_ha"] < ref["lumo_ha"]
    assert ref["sre_ry"] < 1e-8 and ref["states"] >= len(e)
